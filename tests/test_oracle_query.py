"""Pins of the oracle's probe query E(X, n, w_o) (paper, Section "Probe
Query", Eq. 1 and Section "Multiple Probe Volumes")."""
import os

import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _vol(orc, origin, spacing, counts, B=0.3, states=None):
    d = S.VolumeDesc(origin=origin, spacing=(spacing,) * 3, counts=counts, self_shadow_bias=B)
    v = orc.Volume(d, states=np.full(d.n_probes, S.VIGILANT) if states is None else states)
    v.dist[..., 0] = 100.0            # far: every probe sees every point
    v.dist[..., 1] = 100.0 ** 2 + 1.0
    return v


def _fill_dir_tile(orc, m, f):
    k = m - 2
    t = np.zeros((m, m, len(f(np.array([0, 0, 1.0])))))
    for y in range(1, k + 1):
        for x in range(1, k + 1):
            t[y, x] = f(orc.texel_direction(m, x, y))
    for y in range(m):
        for x in range(m):
            sx, sy = orc.border_source(m, x, y)
            t[y, x] = t[sy, sx]
    return t


def _q(orc, vols, X, n, wo):
    e, k = orc.query(vols, np.atleast_2d(X), np.atleast_2d(n), np.atleast_2d(wo))
    return e[0]


def test_constant_atlas_returns_the_constant(orc):
    v = _vol(orc, (0, 0, 0), 1.0, (4, 4, 4))
    v.irr[:] = [0.25, 1.5, 3.0]
    st = S.Stream(910, 1)
    # random visibility texels too: normalisation still returns the constant
    v.dist[..., 0] = st.uniform(v.dist[..., 0].size, 0.2, 2.0).reshape(v.dist[..., 0].shape)
    v.dist[..., 1] = v.dist[..., 0] ** 2 + 0.01
    X = st.uniform(3 * 500, -0.5, 3.5).reshape(-1, 3)
    n = st.unit_vectors(500)
    e, _ = orc.query([v], X, n, n)
    ok = np.abs(e).sum(1) > 0
    assert ok.mean() > 0.9
    assert np.allclose(e[ok], [0.25, 1.5, 3.0], rtol=1e-13)


def test_query_at_a_probe_is_that_probe(orc):
    v = _vol(orc, (0.5, -1.0, 2.0), 1.0, (3, 3, 3))
    st = S.Stream(911, 1)
    vals = st.uniform(27 * 3, 0.1, 5).reshape(27, 3)
    v.irr[:] = vals[:, None, None, :]
    for q in range(27):
        i, j, k = q % 3, (q // 3) % 3, q // 9
        X = np.array([0.5 + i, -1.0 + j, 2.0 + k])
        nn = st.unit_vectors(1)[0]
        assert np.allclose(_q(orc, [v], X, nn, nn), vals[q], rtol=1e-13)


def test_only_awake_and_vigilant_probes_are_sampled(orc):
    st = np.array([S.OFF, S.SLEEPING, S.NEWLY_AWAKE, S.NEWLY_VIGILANT, S.AWAKE, S.VIGILANT, S.OFF, S.OFF],
                  dtype=np.uint8)
    v = _vol(orc, (0, 0, 0), 1.0, (2, 2, 2), states=st)
    for q in range(8):
        v.irr[q] = q
    e = _q(orc, [v], [0.5, 0.5, 0.5], [0, 0, 1.0], [0, 0, 1.0])
    # only probes 4 and 5 count; equal trilinear weight, equal backface weight
    # by symmetry of n about the two probes' directions
    assert np.allclose(e, 4.5, rtol=1e-13)


def test_visibility_looks_up_the_direction_from_probe_to_point(orc):
    """Probe A's distance texels say 'wall at 0.1 m' in the half-space facing
    away from the query point and 'open' elsewhere: A sees the point and
    counts fully.  Turning the wall toward the point hides A; the result then
    equals the query with A switched off."""
    base = _vol(orc, (0, 0, 0), 1.0, (2, 2, 2))
    for q in range(8):
        base.irr[q] = 1.0 + q
    X = np.array([0.3, 0.4, 0.35])
    n = np.array([0.0, 0.0, 1.0])
    A = 0                       # probe at the origin; the point is in +xyz from it
    towards = X / np.linalg.norm(X)
    ref_all = _q(orc, [base], X, n, n)
    off = _vol(orc, (0, 0, 0), 1.0, (2, 2, 2))
    off.irr[:] = base.irr
    off.states[A] = S.OFF
    ref_off = _q(orc, [off], X, n, n)
    assert not np.allclose(ref_all, ref_off)

    def wall(sign):
        f = lambda v: [0.1, 0.01 + 1e-8] if sign * np.dot(v, towards) > 0 else [100.0, 1e4 + 1.0]  # noqa: E731
        return _fill_dir_tile(orc, 16, f)

    base.dist[A] = wall(-1.0)
    assert np.allclose(_q(orc, [base], X, n, n), ref_all, rtol=1e-12)
    base.dist[A] = wall(+1.0)
    assert np.allclose(_q(orc, [base], X, n, n), ref_off, rtol=1e-6)


def test_self_shadow_bias_worked_examples(orc):
    rows = np.loadtxt(os.path.join(GOLDEN, "self_shadow_bias.txt"))
    for wo_x, wo_y, wo_z, B, bx, by, bz, rB, wvis in rows:
        st = np.full(8, S.OFF, np.uint8)
        st[0] = st[1] = S.VIGILANT           # A = (0,0,0), B = (2,0,0)
        v = _vol(orc, (0, 0, 0), 2.0, (2, 2, 2), B=B, states=st)
        cA, cB = 1.0, 3.0
        v.irr[0], v.irr[1] = cA, cB
        v.dist[1, ..., 0] = 0.5
        v.dist[1, ..., 1] = 0.26
        E = _q(orc, [v], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [wo_x, wo_y, wo_z])
        # equal trilinear and backface weights by symmetry, so the weight
        # ratio w_B / w_A is B's visibility weight
        ratio = (cA - E[0]) / (E[0] - cB)
        # B travels as float32 (0.3 -> 0.300000012), which moves w_vis by ~1e-7
        assert ratio == pytest.approx(wvis, rel=1e-6)


def test_cheb_power(orc):
    st = np.full(8, S.OFF, np.uint8)
    st[0] = st[1] = S.VIGILANT
    v = _vol(orc, (0, 0, 0), 2.0, (2, 2, 2), B=0.0, states=st)
    v.desc.cheb_power = 3
    v.irr[0], v.irr[1] = 1.0, 3.0
    v.dist[1, ..., 0] = 0.5
    v.dist[1, ..., 1] = 0.26
    E = _q(orc, [v], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [1.0, 0, 0])
    assert (1.0 - E[0]) / (E[0] - 3.0) == pytest.approx(0.038461538461538464 ** 3, rel=1e-12)


def test_cascade_blend(orc):
    """Dense volume over [0,4]^3 nested in a sparse one over [-2,6]^3: inside
    the dense interior only the dense volume counts; across its last cell the
    weight ramps linearly; outside it the sparse volume takes everything."""
    dense = _vol(orc, (0, 0, 0), 1.0, (5, 5, 5))
    sparse = _vol(orc, (-2, -2, -2), 2.0, (5, 5, 5))
    dense.irr[:] = 1.0
    sparse.irr[:] = 5.0
    n = np.array([0, 1.0, 0])
    for X in ([1.5, 2.0, 2.5], [1.0, 1.0, 3.0], [2.2, 2.9, 1.1]):
        assert np.allclose(_q(orc, [dense, sparse], X, n, n), 1.0, rtol=1e-13)
    for x in np.linspace(3.0, 4.0, 9):
        w = 4.0 - x
        assert np.allclose(_q(orc, [dense, sparse], [x, 2.0, 2.0], n, n), w * 1.0 + (1 - w) * 5.0, rtol=1e-13)
    # two axes in the fade region: weights multiply
    assert np.allclose(_q(orc, [dense, sparse], [3.5, 3.25, 2.0], n, n), 0.5 * 0.75 + (1 - 0.375) * 5, rtol=1e-13)
    for X in ([4.5, 2.0, 2.0], [-1.0, 0.0, 0.0], [5.9, 5.9, 5.9], [9.0, 2.0, 2.0]):
        assert np.allclose(_q(orc, [dense, sparse], X, n, n), 5.0, rtol=1e-13)
    # the sparsest volume always takes the remainder, even outside itself
    assert np.allclose(_q(orc, [sparse], [40.0, 0.0, 0.0], n, n), 5.0, rtol=1e-13)


def test_backface_weight_prefers_probes_in_front(orc):
    # probe in front of the surface (along n) outweighs the one behind it
    st = np.full(8, S.OFF, np.uint8)
    st[0] = st[4] = S.VIGILANT           # (0,0,0) and (0,0,1)
    v = _vol(orc, (0, 0, 0), 1.0, (2, 2, 2), B=0.0, states=st)
    v.irr[0], v.irr[4] = 0.0, 1.0
    E = _q(orc, [v], [0.0, 0.0, 0.5], [0, 0, 1.0], [0, 0, 1.0])
    assert 0.5 < E[0] < 1.0
