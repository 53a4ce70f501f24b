"""Ragged shapes against the FP64 oracle: two volumes whose ray counts (96
and 32) are not multiples of the 64-lane wave, odd probe counts, and four
lights (the room's sun plus three point lights) -- so trace waves straddle
probe and volume boundaries, each wave's shadow slice mixes lights and
probes, and the per-batch slice map, the shadow origins carried by the tasks
and the light-side point-light segments are all exercised; the state step
runs with the room's dynamic box.  Two update frames (ray records, texels,
states) and the query on both volumes."""
import numpy as np
import pytest

from paper_2009_10796_amd import scenes as S
from tests import gpu_helpers as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _workload():
    w = S.config0()
    w.volumes = [
        S.VolumeDesc(origin=(1.3, 1.1, 1.2), spacing=(2.7, 2.9, 2.6), counts=(3, 2, 3), rays_per_probe=96),
        S.VolumeDesc(origin=(0.7, 0.6, 0.9), spacing=(1.55, 1.7, 1.45), counts=(5, 3, 5), rays_per_probe=32),
    ]
    L = w.lights
    w.lights = S.Lights(L.dir_to_light, L.dir_irradiance,
                        np.array([[4.1, 6.3, 3.7], [1.6, 2.2, 6.4], [6.6, 4.4, 1.9]], np.float32),
                        np.array([[8.0, 6.0, 4.0], [3.0, 5.0, 9.0], [6.0, 6.0, 6.0]], np.float32),
                        np.array([0.1, 0.2, 0.3], np.float32))
    return w


def test_ragged_volumes_and_mixed_lights(torch):
    import oracle
    from paper_2009_10796_amd import irf
    w = _workload()
    ctx = irf.build_workload(w)
    osc = oracle.Scene(w.scene)
    ov = [oracle.Volume(d) for d in w.volumes]
    ctx.classify(w.classify_rotations)
    oracle.classify(osc, ov, w.classify_rotations)
    print(f"[ragged] classification differs on {G.copy_states(ctx, ov, torch)} probes", flush=True)
    verdicts = []
    shadow_rays = 0
    for f in (1, 2):
        vs, rep, rec_o, _ = G.frame(torch, ctx, osc, ov, w.lights, w.frame_rotation(f), f"ragged frame {f}")
        verdicts += vs
        shadow_rays += ctx.frame_stats()["shadow_rays"]
        # the first volume ends mid-wave (17 active probes x 96 rays), the frame
        # in a partial wave
        assert len(ctx.ray_records(0)) % 64 != 0 and len(rec_o) % 64 != 0
        for v in range(len(ctx.volumes)):
            assert len(ctx.ray_records(v)) % w.volumes[v].rays_per_probe == 0
    assert shadow_rays > 0
    verdicts += G.queries(torch, ctx, ov, S.surface_points(w.scene, 6000, 0), "ragged")
    G.check(verdicts)
    ctx.close()
