"""Pins of the oracle's convergence refinements (paper, Sections
"Perception-based exponential encoding" and "Fast Convergence Heuristics"):
irradiance texels stored as the new mean to the power 1/gamma and blended in
that encoding; the query decodes each probe's sample to the power gamma/2,
blends, and squares; per-texel thresholds lower the irradiance hysteresis by
0.15 above a change of 0.25 and to 0 above 0.8 (largest per-channel change in
stored units).  Pinned by closed forms on scenes where every quantity is
uniform (no geometry under a sky, the furnace) and by hand-set atlases."""
import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S

G = 5.0


def _desc(gamma=G, thresholds=False, a=0.875, counts=(3, 2, 2), rays=64, **kw):
    return S.VolumeDesc(origin=(0, 0, 0), spacing=(1, 1, 1), counts=counts, rays_per_probe=rays,
                        hysteresis_irr=a, hysteresis_dist=a, irradiance_gamma=gamma, texel_thresholds=thresholds,
                        **kw)


def _frame(orc, sc, v, sky, f):
    orc.update_frame(sc, S.no_lights(sky=sky), [v], S.rotations(0, 1, start_frame=40 + f)[0], records=False)


def _query_all(orc, v, n=200, seed=1):
    st = S.Stream(960, seed)
    X = st.uniform(3 * n, 0.0, 1.0).reshape(-1, 3) * [2.0, 1.0, 1.0]
    nrm = st.unit_vectors(n)
    return orc.query([v], X, nrm, nrm)[0]


def test_encoded_uniform_sky(orc):
    """Converge frame under a uniform sky: every irradiance texel is
    L^(1/gamma); the query decodes to L exactly; distances are unaffected."""
    sc = orc.Scene(S.empty_scene())
    L = np.float32([0.4, 0.9, 1.3]).astype(np.float64)
    v = orc.Volume(_desc())
    _frame(orc, sc, v, L, 0)
    assert np.allclose(v.irr, L ** (1.0 / G), rtol=1e-13)
    dmax = v.desc.resolved_max_distance()
    assert np.allclose(v.dist[..., 0], dmax, rtol=1e-13)
    assert np.allclose(_query_all(orc, v), L, rtol=1e-12)


def _light_to_dark(orc, gamma):
    """Sky L1 for the converge frame, then L0: the stored value follows
    x_k = a x_{k-1} + (1 - a) L0^(1/gamma) and the query returns x_k^gamma."""
    sc = orc.Scene(S.empty_scene())
    L1, L0 = 1.0, 0.01
    a = 0.875
    v = orc.Volume(_desc(gamma=gamma, a=a))
    _frame(orc, sc, v, (L1,) * 3, 0)
    x = L1 ** (1.0 / gamma)
    out = []
    for f in range(1, 12):
        _frame(orc, sc, v, (np.float32(L0),) * 3, f)
        x = a * x + (1 - a) * float(np.float32(L0)) ** (1.0 / gamma)
        assert np.allclose(v.irr, x, rtol=1e-12), f
        E = _query_all(orc, v, n=50, seed=f)
        assert np.allclose(E, x ** gamma, rtol=1e-11), f
        out.append(x ** gamma)
    return out


@pytest.mark.parametrize("gamma", [1.0, G])
def test_light_to_dark_transition_closed_form(orc, gamma):
    _light_to_dark(orc, gamma)


def test_encoding_converges_faster_light_to_dark(orc):
    lin = _light_to_dark(orc, 1.0)
    enc = _light_to_dark(orc, G)
    # every frame after the drop is darker (closer to L0) with the encoding
    assert all(e < l for e, l in zip(enc, lin))
    assert enc[4] < 0.5 * lin[4]


def test_furnace_with_encoding(orc):
    """Closed sphere of emission Le and albedo rho: with the encoding the
    stored value follows x_1 = Le^(1/g), x_k = a x + (1 - a)(Le + rho x^g)^(1/g)
    (a uniform encoded atlas queries to x^g)."""
    Le = np.array([1.0, 2.0, 0.5])
    rho = 0.6
    a = 0.75
    sc = orc.Scene(S.sphere_scene(4.0, 2, emission=Le.tolist(), albedo=rho))
    v = orc.Volume(S.VolumeDesc(origin=(-1, -1, -1), spacing=(1, 1, 1), counts=(3, 3, 3), rays_per_probe=64,
                                hysteresis_irr=a, hysteresis_dist=a, max_distance=20.0, irradiance_gamma=G))
    x = np.zeros(3)
    for f in range(6):
        orc.update_frame(sc, S.no_lights(), [v], S.rotations(0, 1, start_frame=20 + f)[0], records=False)
        x = Le ** (1 / G) if f == 0 else a * x + (1 - a) * (Le + rho * x ** G) ** (1 / G)
        assert np.allclose(v.irr, x, rtol=1e-12), f


def _uniform_blend(orc, old, L, a, gamma, thresholds, d_old=1.0, d_new=3.0):
    """One probe's blend under rays that all carry radiance L and distance
    d_new, from texels old (irradiance) and d_old (mean distance)."""
    n = 64
    omega = orc.sf_directions(n, np.eye(3, dtype=np.float32))
    rgb = np.tile(np.asarray(L, np.float64), (n, 1))
    d = np.full(n, d_new)
    irr = np.zeros((8, 8, 3))
    irr[:] = old
    dist = np.zeros((16, 16, 2))
    dist[..., 0] = d_old
    dist[..., 1] = d_old ** 2
    orc.blend_probe_ex(omega, rgb, d, 50.0, a, a, gamma, thresholds, irr, dist)
    return irr, dist


@pytest.mark.parametrize("change,expect_a", [(0.2, 0.875), (0.5, 0.725), (0.9, 0.0)])
def test_texel_thresholds_levels(orc, change, expect_a):
    old = np.array([0.3, 0.3, 0.3])
    L = old + [0.0, change, 0.0]          # the largest per-channel change decides for all channels
    irr, dist = _uniform_blend(orc, old, L, 0.875, 1.0, True)
    assert np.allclose(irr[1:7, 1:7], expect_a * old + (1 - expect_a) * L, rtol=1e-14)
    # distance texels keep the base hysteresis whatever the change
    assert np.allclose(dist[1:15, 1:15, 0], 0.875 * 1.0 + 0.125 * 3.0, rtol=1e-14)
    # off: the base hysteresis
    irr0, _ = _uniform_blend(orc, old, L, 0.875, 1.0, False)
    assert np.allclose(irr0[1:7, 1:7], 0.875 * old + 0.125 * L, rtol=1e-14)


def test_texel_threshold_floor_and_sign(orc):
    # a small base hysteresis does not go below 0; a drop counts like a rise
    old = np.array([0.9, 0.9, 0.9])
    irr, _ = _uniform_blend(orc, old, old - [0.5, 0.0, 0.0], 0.1, 1.0, True)
    assert np.allclose(irr[1:7, 1:7], old - [0.5, 0.0, 0.0], rtol=1e-14)


def test_texel_thresholds_measure_encoded_change(orc):
    """With the encoding the change is measured in stored units: a linear
    change of 0.19 is an encoded change of 0.327 (> 0.25)."""
    L_old, L_new = 0.01, 0.2
    e_old, e_new = L_old ** (1 / G), L_new ** (1 / G)
    assert L_new - L_old < 0.25 < e_new - e_old < 0.8
    irr, _ = _uniform_blend(orc, np.full(3, e_old), np.full(3, L_new), 0.875, G, True)
    assert np.allclose(irr[1:7, 1:7], 0.725 * e_old + 0.275 * e_new, rtol=1e-13)
    irr, _ = _uniform_blend(orc, np.full(3, e_old), np.full(3, L_new), 0.875, G, False)
    assert np.allclose(irr[1:7, 1:7], 0.875 * e_old + 0.125 * e_new, rtol=1e-13)


def test_query_blends_on_a_gamma_two_curve(orc):
    """Midpoint of a cage edge with the normal across the edge: the two
    probes get equal weights, so E = ((e1^(g/2) + e2^(g/2)) / 2)^2 -- neither
    the linear mean of the decoded values nor the decoded mean."""
    v = orc.Volume(_desc(counts=(2, 2, 2)), states=np.full(8, S.VIGILANT))
    v.dist[..., 0] = 100.0
    v.dist[..., 1] = 100.0 ** 2 + 1.0
    e1, e2 = 0.5, 0.9
    v.irr[:] = 0.0
    v.irr[0] = e1          # probe (0,0,0)
    v.irr[1] = e2          # probe (1,0,0)
    X = np.array([[0.5, 0.0, 0.0]])
    n = np.array([[0.0, 0.0, -1.0]])    # perpendicular to the edge, facing away from the z = 1 probes
    E = orc.query([v], X, n, n)[0][0]
    expect = ((e1 ** 2.5 + e2 ** 2.5) / 2) ** 2
    assert np.allclose(E, expect, rtol=1e-12)
    assert not np.isclose(expect, (e1 ** 5 + e2 ** 5) / 2, rtol=1e-3)
    assert not np.isclose(expect, ((e1 + e2) / 2) ** 5, rtol=1e-3)


def test_threshold_ambiguity_enters_the_sensitivity(orc):
    """A texel whose change sits within float32 rounding of a threshold
    carries the jump between the two outcomes in its sensitivity."""
    sc = orc.Scene(S.empty_scene())
    a = 0.875
    v = orc.Volume(_desc(gamma=1.0, thresholds=True, a=a))
    _frame(orc, sc, v, (0.5, 0.5, 0.5), 0)
    k0 = v.irr_kappa.max()
    # change of exactly 0.25 (+ float32 rounding of the sky)
    _frame(orc, sc, v, (0.75, 0.5, 0.5), 1)
    jump = 0.15 * 0.25
    assert v.irr_kappa.max() * 8 * 2.0 ** -24 >= 0.9 * jump
    # far from a threshold: no jump term
    v2 = orc.Volume(_desc(gamma=1.0, thresholds=True, a=a))
    _frame(orc, sc, v2, (0.5, 0.5, 0.5), 0)
    _frame(orc, sc, v2, (0.6, 0.5, 0.5), 1)
    assert v2.irr_kappa.max() * 8 * 2.0 ** -24 < 1e-5
    assert k0 < 1e3
