"""Pins of the oracle's tracking window and camera-aware volume blending
(paper, Sections "Tracking Windows" and "Multiple Probe Volumes").

The window moves in whole cells when the camera is more than one spacing
from its centre along an axis; surviving probes keep their data at the same
world positions (circular buffer: only the storage phase changes); the
planes that enter are reset and classified; a tracking volume's blend weight
is the per-axis ramp tightened by one cell and centred on the camera, so a
leapfrog does not change what any shaded point sees."""
import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S

ROT = S.rotations(0, 5, start_frame=1000)


def _vol(orc, counts=(5, 3, 4), spacing=1.0, origin=(0.0, 0.0, 0.0), tracking=True):
    d = S.VolumeDesc(origin=origin, spacing=(spacing,) * 3, counts=counts, rays_per_probe=64, tracking=tracking)
    v = orc.Volume(d, states=np.full(d.n_probes, S.VIGILANT))
    v.dist[..., 0] = 100.0            # far: every probe sees every point
    v.dist[..., 1] = 100.0 ** 2 + 1.0
    return v


def _world(v):
    """World position of every storage slot, from the volume's own state."""
    n = np.asarray(v.desc.counts)
    q = np.arange(v.desc.n_probes)
    s = np.stack([q % n[0], (q // n[0]) % n[1], q // (n[0] * n[1])], 1)
    g = (s - v.phase) % n
    return v.origin.astype(np.float64) + g * np.asarray(v.desc.spacing)


def _query(orc, vols, X, n=(0.0, 1.0, 0.0)):
    X = np.atleast_2d(np.asarray(X, np.float64))
    N = np.tile(np.asarray(n, np.float64), (len(X), 1))
    return orc.query(vols, X, N, N)[0]


def test_shift_keeps_surviving_probes_at_their_world_positions(orc):
    sc = orc.Scene(S.empty_scene())
    v = _vol(orc)
    st = S.Stream(970, 1)
    vals = st.uniform(v.desc.n_probes * 3, 0.1, 5.0).reshape(-1, 3)
    v.irr[:] = vals[:, None, None, :]
    before = {tuple(np.round(p, 9)): vals[q] for q, p in enumerate(_world(v))}
    center = np.array([2.0, 1.0, 1.5])
    assert np.allclose(v.camera, center)
    shift = orc.track_volume(sc, v, center + [1.5, -0.2, 0.99], ROT)
    assert list(shift) == [1, 0, 0]
    assert np.allclose(v.origin, [1.0, 0.0, 0.0])
    after = _world(v)
    kept = 0
    for q, p in enumerate(after):
        key = tuple(np.round(p, 9))
        if key in before:
            kept += 1
            assert np.array_equal(v.irr[q, 3, 3], vals[q])          # the slot did not move
            assert np.array_equal(v.irr[q, 3, 3], before[key])      # same probe, same place
            assert v.states[q] == S.VIGILANT
        else:
            # the plane that entered in front: reset and classified (empty space)
            assert p[0] == 1.0 + 4.0
            assert np.all(v.irr[q] == 0.0) and np.all(v.dist[q] == 0.0)
            assert v.states[q] == S.SLEEPING
    assert kept == 4 * 3 * 4
    # queries at surviving probes return their values (the cage follows the phase)
    for q, p in enumerate(after):
        if p[0] < 5.0:
            assert np.allclose(_query(orc, [v], p)[0], vals[q], rtol=1e-13)


def test_negative_shift_and_teleport(orc):
    sc = orc.Scene(S.empty_scene())
    v = _vol(orc)
    v.irr[:] = 1.0
    shift = orc.track_volume(sc, v, [2.0 - 2.5, 1.0, 1.5 + 1.01], ROT)
    assert list(shift) == [-2, 0, 1]
    assert np.allclose(v.origin, [-2.0, 0.0, 1.0])
    assert list(v.phase) == [3, 0, 1]
    w = _world(v)
    fresh = (w[:, 0] < 0.0) | (w[:, 2] > 3.0)
    assert np.all(v.irr[fresh] == 0.0) and np.all(v.irr[~fresh] == 1.0)
    # a jump beyond the window resets every probe
    shift = orc.track_volume(sc, v, [40.0, 1.0, 2.5], ROT)
    assert shift[0] >= 5
    assert np.all(v.irr == 0.0) and np.all(v.states == S.SLEEPING)
    assert abs(v.origin[0] + 2.0 - 40.0) <= 1.0 + 1e-6


def test_new_planes_go_through_the_state_machine(orc):
    # a wall just beyond the window's +x face: the entering plane sees it
    mb = S.MeshBuilder()
    mb.grid_quad((5.6, -1.0, -1.0), (0.0, 0.0, 6.0), (0.0, 4.0, 0.0), 1, 1, material=0)
    sc = orc.Scene(mb.build([[0.5, 0.5, 0.5]], [[0, 0, 0]]))
    v = _vol(orc)
    orc.track_volume(sc, v, [3.5, 1.0, 1.5], ROT)
    w = _world(v)
    front = w[:, 0] == 5.0
    assert np.all(v.states[front] == S.NEWLY_VIGILANT)      # a front face within one spacing
    assert np.all(v.states[~front] == S.VIGILANT)


def test_camera_centred_blend_weight(orc):
    """Dense tracking volume of constant A inside a sparse volume of constant
    B: E = w A + (1 - w) B with w = prod_a clamp(h - |X_a - cam_a| / s, 0, 1),
    h = (n - 1) / 2 - 1."""
    A, B = 2.0, 0.5
    dense = _vol(orc, counts=(7, 7, 7), origin=(0.0, 0.0, 0.0))
    dense.irr[:] = A
    sparse = _vol(orc, counts=(4, 4, 4), spacing=4.0, origin=(-4.0, -4.0, -4.0), tracking=False)
    sparse.irr[:] = B
    c = np.array([3.0, 3.0, 3.0])
    for dx, w in [(1.0, 1.0), (1.5, 0.5), (1.75, 0.25), (2.5, 0.0)]:   # float32-exact points
        E = _query(orc, [dense, sparse], c + [dx, 0.0, 0.0])[0]
        assert np.allclose(E, w * A + (1 - w) * B, rtol=1e-12), dx
    # two axes multiply
    E = _query(orc, [dense, sparse], c + [1.5, -1.75, 0.0])[0]
    assert np.allclose(E, 0.5 * 0.25 * A + (1 - 0.125) * B, rtol=1e-12)
    # the camera moves within its cell: the ramp moves with it (no shift yet)
    sc = orc.Scene(S.empty_scene())
    assert list(orc.track_volume(sc, dense, c + [0.375, 0.0, 0.0], ROT)) == [0, 0, 0]
    E = _query(orc, [dense, sparse], c + [1.5, 0.0, 0.0])[0]
    assert np.allclose(E, 0.875 * A + 0.125 * B, rtol=1e-12)
    # the same point in a non-tracking volume of the same grid: full weight
    static = _vol(orc, counts=(7, 7, 7), origin=(0.0, 0.0, 0.0), tracking=False)
    static.irr[:] = A
    assert np.allclose(_query(orc, [static, sparse], c + [1.5, 0.0, 0.0])[0], A, rtol=1e-12)


def test_leapfrog_does_not_pop(orc):
    """Across a window shift the shaded points see the same probes with
    continuously varying weight: only planes outside the tightened region
    are reinitialised."""
    sc = orc.Scene(S.empty_scene())
    dense = _vol(orc, counts=(7, 7, 7))
    dense.irr[:] = (1.0 + 0.3 * _world(dense)[:, 0])[:, None, None, None]   # varies along x
    sparse = _vol(orc, counts=(4, 4, 4), spacing=4.0, origin=(-4.0, -4.0, -4.0), tracking=False)
    sparse.irr[:] = 0.5
    st = S.Stream(971, 2)
    X = st.uniform(3 * 400, 0.0, 7.0).reshape(-1, 3)
    c = np.array([3.0, 3.0, 3.0])
    orc.track_volume(sc, dense, c + [0.999, 0.0, 0.0], ROT)
    E1 = _query(orc, [dense, sparse], X)
    assert list(orc.track_volume(sc, dense, c + [1.001, 0.0, 0.0], ROT)) == [1, 0, 0]
    E2 = _query(orc, [dense, sparse], X)
    # the weights moved by 0.002 of a cell: E moves by at most that fraction of |A - B|
    assert np.max(np.abs(E2 - E1)) <= 0.002 * (1.0 + 0.3 * 7.0) + 1e-12
