"""The query-stage tolerance of the GPU parity tests is tight enough to see
a texel fetched from the wrong place: on the oracle's own converged room
(atlases rounded to float16, as the half-atlas GPU test stores them), the
two texels of every horizontal pair of a tile row are swapped -- in the
irradiance tiles, then in the distance tiles -- and the oracle's query of
the planted atlas must fall outside the tolerance for many points.  (A
swapped pair is what a wrong wide load of adjacent texels would produce.)"""
import numpy as np

from paper_2009_10796_amd import scenes as S
from tests import parity as P


def _swap_pairs(a):
    s = a.copy()
    s[:, :, 0::2], s[:, :, 1::2] = a[:, :, 1::2].copy(), a[:, :, 0::2].copy()
    return s


def test_swapped_texel_pairs_fail_the_query_tolerance():
    import oracle
    w = S.config0(n_queries=20000)
    for d in w.volumes:
        d.atlas_f16 = True
    osc = oracle.Scene(w.scene)
    ov = [oracle.Volume(d) for d in w.volumes]
    oracle.classify(osc, ov, w.classify_rotations)
    for f in (1, 2):
        oracle.update_frame(osc, w.lights, ov, w.frame_rotation(f), records=False)
    o = ov[0]
    irr = o.irr.astype(np.float16).astype(np.float64)
    dist = o.dist.astype(np.float16).astype(np.float64)

    def query(i, d):
        v = oracle.Volume(w.volumes[0], states=o.states)
        v.irr[:] = i
        v.dist[:] = d
        return oracle.query([v], w.queries.pos, w.queries.nrm, w.queries.view)

    eo, ko = query(irr, dist)
    assert P.compare("unchanged", eo, eo, ko).ok
    for planted in (query(_swap_pairs(irr), dist)[0], query(irr, _swap_pairs(dist))[0]):
        v = P.compare("planted", planted, eo, ko)
        assert v.fail > 0.1 * eo.size, v.line()
