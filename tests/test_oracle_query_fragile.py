"""The oracle's float32 sensitivity of a query whose every weight is
undetermined in float32 (Section "Probe Query": weights normalised by their
sum; zero when no probe carries weight).

One sampled probe of a 2x2x2 volume, queried beyond its distance clamp, so
its weight is the one-sided Chebyshev bound var / (var + (r - mu)^2).  With
the stored mean square at mu^2 (1 + 1e-9) the variance lies below the
float32 resolution of mu2 - mu^2: float32 may find it zero, the weight sum
zero and the query zero, while the exact result is the probe's irradiance
(the normalisation removes the tiny weight).  The oracle's kappa must then
cover the whole value (8 u kappa >= |E|).  With mu^2 (1 + 1e-3) the
variance is resolved and kappa stays a small multiple of |E|."""
import numpy as np

from paper_2009_10796_amd import scenes as S

U32 = 2.0 ** -24


def _query(rel_excess):
    import oracle
    d = S.VolumeDesc(origin=(0.0, 0.0, 0.0), spacing=(1.0, 1.0, 1.0), counts=(2, 2, 2), rays_per_probe=64)
    states = np.zeros(8, np.uint8)
    states[1] = S.VIGILANT                       # the probe at (1, 0, 0)
    v = oracle.Volume(d, states=states)
    mu = d.resolved_max_distance()
    v.irr[1] = np.array([1.0, 2.0, 3.0])
    v.dist[1, ..., 0] = mu
    v.dist[1, ..., 1] = mu * mu * (1.0 + rel_excess)
    X = np.array([[4.0, 0.0, 0.0]], np.float32)   # clamped cage: all weight on the x = 1 plane
    n = np.array([[-1.0, 0.0, 0.0]], np.float32)  # facing the probe
    E, k = oracle.query([v], X, n, n)
    return E[0], k[0]


def test_fragile_only_weight_covers_a_zero_result():
    E, k = _query(1e-9)
    assert np.allclose(E, [1.0, 2.0, 3.0], rtol=1e-9)
    assert np.all(8 * U32 * k >= np.abs(E))


def test_resolved_variance_keeps_kappa_small():
    E, k = _query(1e-3)
    assert np.allclose(E, [1.0, 2.0, 3.0], rtol=1e-9)
    assert np.all(8 * U32 * k < 1e-3 * np.abs(E))
