"""Pins of the oracle's ray directions and nearest-hit search.

Probe rays follow a spherical-Fibonacci pattern with a random rotation per
frame (paper, Section "Probe Update").  The nearest hit is a plain minimum
over triangles; the oracle's own BVH is only an accelerator and is pinned to
brute force here, and brute force is pinned to analytic geometry.
"""
import math

import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S

PHI = (1 + 5 ** 0.5) / 2


def test_sf_closed_form_and_uniformity(orc):
    I = np.eye(3, dtype=np.float32)
    for n in (64, 192, 256, 1024):
        w = orc.sf_directions(n, I)
        i = np.arange(n)
        assert np.allclose(w[:, 2], 1 - (2 * i + 1) / n, atol=1e-15)          # equal-area bands
        assert np.allclose(np.linalg.norm(w, axis=1), 1.0, atol=1e-14)
        assert abs(w[:, 2].sum()) < 1e-11
        # azimuth advances by the golden angle 2*pi*(phi - 1)
        az = np.arctan2(w[:, 1], w[:, 0])
        step = np.mod(np.diff(az), 2 * np.pi)
        assert np.allclose(step, np.mod(2 * np.pi * (PHI - 1), 2 * np.pi), atol=1e-9)
        # quadrature of low-order moments of the uniform sphere
        assert np.allclose(w.mean(0), 0.0, atol=2.0 / n)
        assert abs((w[:, 2] ** 2).mean() - 1 / 3) < 1.0 / n
        assert abs((w[:, 0] ** 2).mean() - 1 / 3) < 4.0 / n


def test_rotation_applies_to_the_pattern(orc):
    R = S.rotations(0, 1)[0]
    I = np.eye(3, dtype=np.float32)
    base = orc.sf_directions(64, I)
    rot = orc.sf_directions(64, R)
    assert np.allclose(rot, base @ R.reshape(3, 3).astype(np.float64).T, atol=1e-14)


def test_room_walls_analytic(orc):
    """Rays from inside the closed 8 m room hit the walls where the slab
    distance says, when nothing else is in the way."""
    mb = S.MeshBuilder()
    mb.box((0, 0, 0), (8, 8, 8), material=0, inward=True)
    sc = orc.Scene(mb.build([[0.5] * 3], [[0, 0, 0]]))
    o = np.array([2.3, 5.1, 3.7])
    dirs = S.Stream(903, 1).unit_vectors(400)
    hits = sc.trace(np.repeat(o[None], len(dirs), 0), dirs)
    t_exp = np.min(np.where(dirs > 0, (8 - o) / np.where(dirs == 0, 1, dirs),
                            np.where(dirs < 0, (0 - o) / np.where(dirs == 0, 1, dirs), np.inf)), axis=1)
    assert np.all(hits["tri"] >= 0)
    assert np.allclose(hits["t"], t_exp, rtol=1e-13)


def test_bvh_equals_brute_force(orc):
    soup = S.random_triangle_soup(600)
    sc = orc.Scene(soup)
    st = S.Stream(904, 1)
    o = st.uniform(3 * 3000, -5, 5).reshape(-1, 3)
    d = st.unit_vectors(3000)
    for static_only in (False, True):
        a = sc.trace(o, d, static_only=static_only)
        b = sc.trace(o, d, static_only=static_only, brute=True)
        assert np.array_equal(a["tri"], b["tri"])
        assert np.array_equal(a["t"], b["t"])
        assert np.array_equal(a["flags"], b["flags"])
        assert (a["tri"] >= 0).mean() > 0.3
    # the static-only trace never returns a dynamic triangle
    a = sc.trace(o, d, static_only=True)
    hit = a["tri"] >= 0
    assert np.all(soup.tri_object[a["tri"][hit]] == 0)


def test_closed_sphere_is_watertight(orc):
    sc = orc.Scene(S.sphere_scene(radius=3.0, subdiv=3))
    st = S.Stream(905, 1)
    o = st.uniform(3 * 2000, -1.5, 1.5).reshape(-1, 3)
    d = st.unit_vectors(2000)
    h = sc.trace(o, d)
    assert np.all(h["tri"] >= 0)
    # the hit point is on the tessellated sphere: between inscribed and circumscribed radii
    X = o + h["t"][:, None] * d
    r = np.linalg.norm(X, axis=1)
    assert np.all(r <= 3.0 + 1e-12) and np.all(r >= 3.0 * 0.98)


def test_flags_mark_edge_hits(orc):
    # two triangles sharing the edge x = 0 of a unit square in the plane z = 0
    verts = np.array([[-1, -1, 0], [0, -1, 0], [0, 1, 0], [-1, 1, 0], [1, -1, 0], [1, 1, 0]], np.float32)
    idx = np.array([[0, 1, 2], [0, 2, 3], [1, 4, 5], [1, 5, 2]], np.uint32)
    sc = orc.Scene(S.Scene(verts, idx, np.zeros(4, np.uint32), np.zeros(4, np.uint32),
                           np.full((1, 3), 0.5, np.float32), np.zeros((1, 3), np.float32)))
    down = np.array([[0, 0, -1.0]])
    # exactly on the shared edge: a hit, flagged as grazing and as a tie
    h = sc.trace(np.array([[0.0, 0.3, 1.0]]), down)[0]
    assert h["tri"] >= 0 and h["flags"] & orc.F_GRAZE and h["flags"] & orc.F_TIE
    assert h["t"] == 1.0
    # well inside one triangle: unflagged
    h = sc.trace(np.array([[0.5, -0.2, 1.0]]), down)[0]
    assert h["flags"] == 0 and h["t"] == 1.0
    # just outside the outer edge: a miss, flagged as a near miss
    h = sc.trace(np.array([[1.0 + 1e-6, 0.0, 1.0]]), down)[0]
    assert h["tri"] < 0 and h["flags"] & orc.F_NEARMISS
    # far outside: a clean miss
    h = sc.trace(np.array([[3.0, 0.0, 1.0]]), down)[0]
    assert h["tri"] < 0 and h["flags"] == 0


def test_nearest_of_stacked_planes(orc):
    # parallel planes at z = 0, 1, 2 (front +z); a ray down from z = 5 hits z = 2 first
    mb = S.MeshBuilder()
    for z in (0.0, 1.0, 2.0):
        mb.grid_quad((-4, -4, z), (8, 0, 0), (0, 8, 0), 3, 3, material=0)
    sc = orc.Scene(mb.build([[0.5] * 3], [[0, 0, 0]]))
    st = S.Stream(906, 1)
    n = 500
    o = np.column_stack([st.uniform(n, -1, 1), st.uniform(n, -1, 1), np.full(n, 5.0)])
    d = np.column_stack([st.uniform(n, -0.3, 0.3), st.uniform(n, -0.3, 0.3), -np.ones(n)])
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    h = sc.trace(o, d)
    assert np.allclose(h["t"], 3.0 / -d[:, 2], rtol=1e-13)
    # from z = 1.5 upward the z = 2 plane is hit from behind
    h = sc.trace(np.array([[0.1, 0.2, 1.5]]), np.array([[0, 0, 1.0]]))[0]
    assert h["t"] == pytest.approx(0.5, abs=1e-15)
