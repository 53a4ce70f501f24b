"""Pins of the oracle's probe relocation (paper, Section "Probe Position
Adjustment").  The geometry of each case is solved here independently
(rays against axis-aligned walls and a single quad, in numpy), and the
optimizer's move is checked by what the section says it does: through the
closest backface to the edge of the allowed offset box, or a bounded step
toward the farthest front face, or no move."""
import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S

SP = 10.0          # spacing: the other probes of the 2x2x2 volume are far away


def _setup(orc, mb, rays=256):
    sc = orc.Scene(mb.build([[0.5, 0.5, 0.5]], [[0, 0, 0]]))
    d = S.VolumeDesc(origin=(0, 0, 0), spacing=(SP, SP, SP), counts=(2, 2, 2), rays_per_probe=rays)
    return sc, orc.Volume(d)


def _rays(orc, n, R):
    return orc.sf_directions(n, R)


def _box_exit(w, lo, hi, p=np.zeros(3)):
    """Distance from p (inside the box) to the box boundary along each ray."""
    t = np.full(len(w), np.inf)
    for a in range(3):
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = np.where(w[:, a] > 0, (hi[a] - p[a]) / w[:, a], np.where(w[:, a] < 0, (lo[a] - p[a]) / w[:, a], np.inf))
        t = np.minimum(t, ta)
    return t


R0 = S.rotations(0, 5, start_frame=1010)


def test_probe_inside_a_box_moves_through_the_closest_backface(orc):
    lo, hi = np.array([-0.3, -1.0, -1.0]), np.array([1.0, 1.0, 1.0])
    mb = S.MeshBuilder()
    mb.box(lo, hi, material=0)               # outward faces: all backfaces from inside
    sc, v = _setup(orc, mb)
    limit = 0.05                               # 0.5 m per axis
    amb = orc.optimize_offsets(sc, v, R0[:1], offset_limit=limit)
    assert amb[0] == 0
    w = _rays(orc, 256, R0[0])
    t = _box_exit(w, lo, hi)
    r = int(np.argmin(t))
    off = v.offsets[0].astype(np.float64)
    # along the ray to the closest backface ...
    assert np.allclose(off / np.linalg.norm(off), w[r], atol=1e-6)
    # ... past the backface (outside the box) ...
    assert np.linalg.norm(off) > t[r]
    assert np.any(off < lo) or np.any(off > hi)
    # ... to the edge of the offset box, less 1e-3 of the scale
    lim = limit * SP
    s = np.linalg.norm(off) / t[r]
    assert np.isclose(np.max(np.abs(off)) + 1e-3 * np.max(np.abs(w[r] * t[r])), lim, rtol=1e-6)
    assert s > 1


def test_probe_that_cannot_get_through_stays(orc):
    lo, hi = np.array([-0.6, -1.0, -1.0]), np.array([1.0, 1.0, 1.0])
    mb = S.MeshBuilder()
    mb.box(lo, hi, material=0)
    sc, v = _setup(orc, mb)
    orc.optimize_offsets(sc, v, R0[:1], offset_limit=0.05)   # 0.5 m < 0.6 m to the nearest wall
    assert np.all(v.offsets[0] == 0.0)


def _quad_hits(w, o, u, vv, p=np.zeros(3)):
    """Front-face hits of rays from p on the parallelogram o + a u + b v
    (front side u x v); inf where missed or seen from behind."""
    n = np.cross(u, vv)
    den = w @ n
    with np.errstate(divide="ignore", invalid="ignore"):
        t = ((o - p) @ n) / den
    X = p + t[:, None] * w
    M = np.stack([u, vv], 1)
    ab = np.linalg.lstsq(M, (X - o).T, rcond=None)[0].T
    ok = (den < 0) & (t > 0) & (ab[:, 0] >= 0) & (ab[:, 0] <= 1) & (ab[:, 1] >= 0) & (ab[:, 1] <= 1)
    return np.where(ok, t, np.inf)


def test_probe_near_a_wall_steps_toward_the_farthest_front_face(orc):
    # a 3 x 3 m wall 0.3 m in front of the probe, facing it (+x side)
    o, u, vv = np.array([0.3, -1.5, -1.5]), np.array([0.0, 0.0, 3.0]), np.array([0.0, 3.0, 0.0])
    assert np.cross(u, vv)[0] < 0     # front side faces the probe at the origin
    mb = S.MeshBuilder()
    mb.grid_quad(o, u, vv, 1, 1, material=0)
    sc, v = _setup(orc, mb)
    amb = orc.optimize_offsets(sc, v, R0[:1], offset_limit=0.45)
    assert amb[0] == 0
    w = _rays(orc, 256, R0[0])
    t = _quad_hits(w, o, u, vv)
    hit = np.isfinite(t)
    rf = int(np.argmax(np.where(hit, t, -1)))
    rc = int(np.argmin(t))
    assert np.dot(w[rf], w[rc]) <= 0.5          # the wall spans more than 60 degrees
    expect = min(0.2, t[rf]) * w[rf]
    assert np.allclose(v.offsets[0], expect, atol=1e-6)


def test_probe_seeing_one_small_surface_stays(orc):
    # a 0.4 m square 3 m away: every hit within a narrow cone
    o, u, vv = np.array([3.0, -0.2, -0.2]), np.array([0.0, 0.0, 0.4]), np.array([0.0, 0.4, 0.0])
    mb = S.MeshBuilder()
    mb.grid_quad(o, u, vv, 1, 1, material=0)
    sc, v = _setup(orc, mb, rays=1024)
    w = _rays(orc, 1024, R0[0])
    t = _quad_hits(w, o, u, vv)
    assert np.isfinite(t).sum() >= 2
    orc.optimize_offsets(sc, v, R0[:1], offset_limit=0.45)
    assert np.all(v.offsets[0] == 0.0)


def test_empty_scene_and_dynamic_geometry_do_not_move_probes(orc):
    sce = orc.Scene(S.empty_scene())
    v = orc.Volume(S.VolumeDesc(origin=(0, 0, 0), spacing=(1, 1, 1), counts=(2, 2, 2), rays_per_probe=64))
    amb = orc.optimize_offsets(sce, v, R0, offset_limit=0.45)
    assert np.all(v.offsets == 0.0) and np.all(amb == 0)
    # a box that is a dynamic object: not seen by the optimizer
    mb = S.MeshBuilder()
    mb.box((-0.3, -1, -1), (1, 1, 1), material=0, obj=1)
    sc, v = _setup(orc, mb)
    orc.optimize_offsets(sc, v, R0[:1], offset_limit=0.05)
    assert np.all(v.offsets == 0.0)


def test_five_iterations_leave_the_probe_outside_and_in_bounds(orc):
    lo, hi = np.array([-0.3, -1.0, -1.0]), np.array([1.0, 1.0, 1.0])
    mb = S.MeshBuilder()
    mb.box(lo, hi, material=0)
    sc, v = _setup(orc, mb)
    orc.optimize_offsets(sc, v, R0, offset_limit=0.05)
    off = v.offsets[0].astype(np.float64)
    assert np.any(off < lo) or np.any(off > hi)
    assert np.all(np.abs(v.offsets) <= 0.05 * SP + 1e-6)


def test_relocation_reduces_off_probes_in_the_city(orc):
    """City volume: probes inside buildings see backfaces and are classified
    Off; relocation moves those within reach of a wall out."""
    w = S.config1(gbuffer=False)
    sc = orc.Scene(w.scene)
    before = orc.Volume(w.volumes[0])
    orc.classify(sc, [before], w.classify_rotations)
    after = orc.Volume(w.volumes[0])
    amb = orc.optimize_offsets(sc, after, S.rotations(1, 5, start_frame=1010), offset_limit=0.45)
    orc.classify(sc, [after], w.classify_rotations)
    n_off_before = int((before.states == S.OFF).sum())
    n_off_after = int((after.states == S.OFF).sum())
    print(f"Off probes: {n_off_before} -> {n_off_after}; ambiguous {int((amb != 0).sum())}")
    assert n_off_after < n_off_before
    assert np.all(np.abs(after.offsets) <= 0.45 + 1e-6)
