"""Pins of the oracle's octahedral map, texel layout and tile sampling.

The probes store spherical functions in octahedral tiles (Cigolle et al.
2014), 8x8 irradiance and 16x16 distance with a one-texel border for
bilinear filtering (paper, Table 2 and Section "Probe Update Shader
Optimization").  These tests check the oracle against closed forms of the
map and against the geometry of the octahedral seam, not against itself.
"""
import numpy as np
import pytest

from paper_2009_10796_amd.scenes import Stream


def _rand_dirs(n, seed=7):
    return Stream(900, seed).unit_vectors(n)


def test_encode_decode_round_trip(orc):
    dirs = list(_rand_dirs(500)) + [np.array(v, float) for v in
                                     [(1, 0, 0), (0, 1, 0), (0, 0, 1), (0, 0, -1), (-1, 0, 0), (0, -1, 0),
                                      (1, 1, 0), (1, -1, -1e-12), (0.3, -0.2, -0.9)]]
    for v in dirs:
        v = v / np.linalg.norm(v)
        p = orc.oct_encode(v)
        assert np.all(np.abs(p) <= 1.0)
        assert np.allclose(orc.oct_decode(p), v, atol=1e-14)


def test_upper_hemisphere_is_the_inner_diamond(orc):
    # closed form: for z >= 0 the map is the L1-normalised (x, y)
    for v in _rand_dirs(200, 8):
        v[2] = abs(v[2])
        p = orc.oct_encode(v)
        l1 = np.abs(v).sum()
        assert np.allclose(p, v[:2] / l1, atol=1e-15)
        assert abs(p).sum() <= 1 + 1e-15


def test_seam_fold_identities(orc):
    # the square's edges fold onto themselves: (a, +-1) ~ (-a, +-1), (+-1, b) ~ (+-1, -b)
    for a in np.linspace(-1, 1, 17):
        for s in (-1.0, 1.0):
            assert np.allclose(orc.oct_decode([a, s]), orc.oct_decode([-a, s]), atol=1e-15)
            assert np.allclose(orc.oct_decode([s, a]), orc.oct_decode([s, -a]), atol=1e-15)
    # all four corners are the south pole
    for c in [(-1, -1), (-1, 1), (1, -1), (1, 1)]:
        assert np.allclose(orc.oct_decode(c), [0, 0, -1], atol=1e-15)


def _wrap(p):
    """Continuation of the octahedral square across its seam: leaving through
    the edge y = +-1 re-enters mirrored in x; leaving through x = +-1 re-enters
    mirrored in y.  Derived from the fold identities above."""
    x, y = p
    if y > 1:
        x, y = -x, 2 - y
    elif y < -1:
        x, y = -x, -2 - y
    if x > 1:
        x, y = 2 - x, -y
    elif x < -1:
        x, y = -2 - x, -y
    return x, y


@pytest.mark.parametrize("m", [8, 16])
def test_border_cells_hold_the_cell_across_the_seam(orc, m):
    k = m - 2
    centre = lambda c: 2.0 * ((c - 1) + 0.5) / k - 1.0  # noqa: E731  (cell index -> square coordinate)
    for y in range(m):
        for x in range(m):
            sx, sy = orc.border_source(m, x, y)
            if 1 <= x <= k and 1 <= y <= k:
                assert (sx, sy) == (x, y)
                continue
            assert 1 <= sx <= k and 1 <= sy <= k
            wx, wy = _wrap((centre(x), centre(y)))
            assert np.isclose(wx, centre(sx), atol=1e-12) and np.isclose(wy, centre(sy), atol=1e-12), (x, y)


@pytest.mark.parametrize("m", [8, 16])
def test_texel_directions_are_decoded_cell_centres(orc, m):
    k = m - 2
    seen = []
    for y in range(1, k + 1):
        for x in range(1, k + 1):
            v = orc.texel_direction(m, x, y)
            assert np.isclose(np.linalg.norm(v), 1.0, atol=1e-15)
            p = orc.oct_encode(v)
            assert np.allclose(p, [2 * (x - 0.5) / k - 1, 2 * (y - 0.5) / k - 1], atol=1e-14)
            seen.append(v)
    # the interior covers the sphere symmetrically
    assert np.allclose(np.mean(seen, axis=0), 0.0, atol=1e-12)


def _filled_tile(orc, m, f):
    k = m - 2
    tile = np.zeros((m, m, 1))
    for y in range(1, k + 1):
        for x in range(1, k + 1):
            tile[y, x, 0] = f(orc.texel_direction(m, x, y))
    for y in range(m):
        for x in range(m):
            sx, sy = orc.border_source(m, x, y)
            tile[y, x, 0] = tile[sy, sx, 0]
    return tile


@pytest.mark.parametrize("m", [8, 16])
def test_sampling_a_texel_centre_returns_the_texel(orc, m):
    k = m - 2
    tile = _filled_tile(orc, m, lambda v: 0)
    tile[..., 0] = Stream(901, m).uniform(m * m).reshape(m, m)
    for y in range(1, k + 1):
        for x in range(1, k + 1):
            assert orc.sample_tile(tile, orc.texel_direction(m, x, y))[0] == pytest.approx(tile[y, x, 0], abs=1e-12)


@pytest.mark.parametrize("m", [8, 16])
def test_bilinear_is_continuous_across_the_seam(orc, m):
    """With the border filled by the seam rule, the interpolated field is
    continuous on the sphere: two directions just either side of a seam give
    the same sample in the limit.  A border that is not the mirrored cell
    (for example clamp-to-edge) leaves a jump of the size of the data."""
    tile = _filled_tile(orc, m, lambda v: 0)
    tile[..., 0] = Stream(902, m).uniform(m * m).reshape(m, m)
    for y in range(m):
        for x in range(m):
            sx, sy = orc.border_source(m, x, y)
            tile[y, x, 0] = tile[sy, sx, 0]
    d = 1e-9
    for a in np.linspace(-0.97, 0.97, 23):
        for s in (-1.0, 1.0):
            # across the edge y = s: (a, s - s d) and (-a, s - s d)
            v1 = orc.oct_decode([a, s * (1 - d)])
            v2 = orc.oct_decode([-a, s * (1 - d)])
            assert np.linalg.norm(v1 - v2) < 1e-6
            assert abs(orc.sample_tile(tile, v1)[0] - orc.sample_tile(tile, v2)[0]) < 1e-6
            # across the edge x = s
            v1 = orc.oct_decode([s * (1 - d), a])
            v2 = orc.oct_decode([s * (1 - d), -a])
            assert abs(orc.sample_tile(tile, v1)[0] - orc.sample_tile(tile, v2)[0]) < 1e-6
    # near the south pole all four corners meet
    vals = [orc.sample_tile(tile, orc.oct_decode([sx * (1 - d), sy * (1 - d)]))[0]
            for sx in (-1, 1) for sy in (-1, 1)]
    assert max(vals) - min(vals) < 1e-6


def test_sampling_clamps_inside_the_tile(orc):
    # every tap stays inside [0, m-1]: sampling a tile whose border is NaN-free
    # and whose interior is constant returns the constant everywhere
    for m in (8, 16):
        tile = np.full((m, m, 2), 3.25)
        for v in list(_rand_dirs(300, 10)) + [np.array([0, 0, -1.0]), np.array([1.0, 0, 0])]:
            assert np.allclose(orc.sample_tile(tile, v), 3.25, atol=1e-14)
