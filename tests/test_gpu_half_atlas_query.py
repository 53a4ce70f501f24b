"""Query stage on half-precision atlases against the FP64 oracle.

The oracle converges the probes (classification, two update frames); its
atlases, rounded to float16, are stored in the GPU's half atlases and given
back to a fresh oracle volume as the same rounded values, so both sides
query identical texels.  The GPU then reads each bilinear texel pair of a
tile row with one wide load (a half4 irradiance pair as 16 bytes, a half2
distance pair as 8), which the float32-atlas tests do not reach.  Room
(random points, random normals and views: every texel pair of the tiles)
with linear and with perceptually encoded irradiance, and the full city
G-buffer with linear irradiance.  Tolerance as in the float32 query stage."""
import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S
from tests import gpu_helpers as G
from tests import parity as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("name,gamma", [("room", 1.0), ("room", 5.0), ("city", 1.0)])
def test_half_atlas_query_stage(torch, name, gamma):
    import oracle
    from paper_2009_10796_amd import irf
    w = S.config0(n_queries=20000) if name == "room" else S.config1()
    for d in w.volumes:
        d.atlas_f16 = True
        d.irradiance_gamma = gamma
    osc = oracle.Scene(w.scene)
    ov = [oracle.Volume(d) for d in w.volumes]
    oracle.classify(osc, ov, w.classify_rotations)
    for f in (1, 2):
        oracle.update_frame(osc, w.lights, ov, w.frame_rotation(f), records=False)
    o = ov[0]
    irr16 = o.irr.astype(np.float16)
    dist16 = o.dist.astype(np.float16)
    assert np.isfinite(irr16).all() and np.isfinite(dist16).all()
    ctx = irf.build_workload(w)
    gv = ctx.volumes[0]
    assert gv.irradiance.dtype == torch.float16 and gv.distance.dtype == torch.float16
    gv.irradiance[..., :3].copy_(torch.from_numpy(irr16))
    gv.distance.copy_(torch.from_numpy(dist16))
    gv.states.copy_(torch.from_numpy(o.states))
    o16 = oracle.Volume(w.volumes[0], states=o.states)
    o16.irr[:] = irr16.astype(np.float64)
    o16.dist[:] = dist16.astype(np.float64)
    q = w.queries
    sampled = np.isin(o.states, [S.AWAKE, S.VIGILANT]).sum()
    print(f"[half atlas] {name} gamma={gamma}: {q.n} queries, {sampled} sampled probes of {len(o.states)}",
          flush=True)
    assert sampled > 0
    e = ctx.query_irradiance(*(torch.from_numpy(a).cuda() for a in (q.pos, q.nrm, q.view))).cpu().numpy()
    eo, ko = oracle.query([o16], q.pos, q.nrm, q.view)
    nz = int((np.abs(eo).max(1) > 0).sum())
    print(f"[half atlas] {name} gamma={gamma}: {nz} of {len(e)} with irradiance", flush=True)
    assert nz > 0.5 * len(e)
    G.check([P.compare(f"half atlas {name} gamma={gamma} query stage", e, eo, ko)])
    ctx.close()
